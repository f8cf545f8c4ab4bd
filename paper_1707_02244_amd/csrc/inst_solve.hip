// Persistent-solver instantiation for one size N = 2^CS_LOGN (complex points,
// n = 2N reals), untraced (CS_TRACE = 0) or with the objective trace
// (CS_TRACE = 1).  Odd log2 N: N2 = 2 N1, two row pairs per workgroup; even:
// N2 = 4 N1, one row pair per workgroup.
#include "launch.hpp"
#include "solve_persistent.hpp"

#ifndef CS_LOGN
#error "compile with -DCS_LOGN=<log2 of the complex length>"
#endif
#ifndef CS_TRACE
#define CS_TRACE 0
#endif

namespace cs {

namespace {
constexpr int kLogN = CS_LOGN;
constexpr int kN1 = (kLogN % 2) ? (1 << ((kLogN - 1) / 2)) : (1 << (kLogN / 2 - 1));
constexpr int kN2 = (1 << kLogN) / kN1;
constexpr int kAI = (kLogN % 2) ? 2 : 1;
constexpr bool kTR = CS_TRACE != 0;

template <int D2, int ALG>
const void* kernel_ptr() {
  if constexpr (kN2 / D2 >= 2) return reinterpret_cast<const void*>(&k_solve<kN1, kN2, D2, kAI, ALG, kTR>);
  else return nullptr;
}

const void* pick(int alg, int d2) {
  switch (d2) {
    case 1: return alg ? kernel_ptr<1, 1>() : kernel_ptr<1, 0>();
    case 2: return alg ? kernel_ptr<2, 1>() : kernel_ptr<2, 0>();
    case 4: return alg ? kernel_ptr<4, 1>() : kernel_ptr<4, 0>();
    case 8: return alg ? kernel_ptr<8, 1>() : kernel_ptr<8, 0>();
    default: return nullptr;
  }
}
}  // namespace

template <>
hipError_t launch_solve<CS_LOGN, kTR>(int alg, int d2, const SolveArgs& a, hipStream_t s) {
  const void* f = pick(alg, d2);
  if (!f) return hipErrorInvalidValue;
  SolveArgs copy = a;
  void* params[] = {&copy};
  return hipLaunchCooperativeKernel(f, dim3(kN2 / kColsPerBlock), dim3(kPThreads), params, 0, s);
}

template <>
int solve_blocks_per_cu<CS_LOGN, kTR>(int alg, int d2) {
  const void* f = pick(alg, d2);
  if (!f) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kPThreads, 0) != hipSuccess) return 0;
  return nb;
}

}  // namespace cs
