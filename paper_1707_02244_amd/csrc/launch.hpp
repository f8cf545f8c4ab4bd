// Host-side launchers for the kernel templates.  Each size is instantiated in
// its own translation unit (inst_passA.hip / inst_passB.hip compiled once per
// length with -DCS_LEN=<L>) so the build parallelises.
#pragma once
#include <hip/hip_runtime.h>
#include "kernels.hpp"

namespace cs {

template <int N2>
hipError_t launch_passA(int op, int d2, int grid, const PassAArgs& a, hipStream_t s);

template <int N1>
hipError_t launch_passB(int mode, int grid, const PassBArgs& a, hipStream_t s);

}  // namespace cs
