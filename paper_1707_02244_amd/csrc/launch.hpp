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

struct CpArgs;
// circulant ADMM with an arbitrary row set (cpadmm.hpp): row pass over row
// pairs, column pass over column blocks (last: write the outputs)
template <int N2>
hipError_t launch_cp_row(int grid, const CpArgs& a, hipStream_t s);
template <int N1>
hipError_t launch_cp_col(int last, int grid, const CpArgs& a, hipStream_t s);

struct UStride;
// batched (grid y = signal) row / column passes for the unrolled solver
template <int N2>
hipError_t launch_urow(int op, int d2, int grid, int batch, const PassAArgs& a, const UStride& st,
                       hipStream_t s);
template <int N1>
hipError_t launch_ucol(int mode, int grid, int batch, const PassBArgs& a, const UStride& st, hipStream_t s);

struct SolveArgs;
// persistent solver for N = 2^LOGN complex points (inst_solve.hip); TR: the
// instance that also writes the objective trace's partial sums
template <int LOGN, bool TR>
hipError_t launch_solve(int alg, int d2, const SolveArgs& a, hipStream_t s);
template <int LOGN, bool TR>
int solve_blocks_per_cu(int alg, int d2);

// persistent batched solver, ALG 0: ISTA, 1: ADMM (inst_bpersist.hip): the
// kernel (launched cooperatively with one PBatchArgs argument) and how many
// of its workgroups fit on one CU
template <int ALG>
const void* batch_persist_kernel();
template <int ALG>
int batch_persist_blocks_per_cu();

struct Col2Args;
struct Row2Args;
// 2-D path: column pass over R-point columns, row pass over H-point rows
// (inst2d_col.hip / inst2d_row.hip)
template <int R>
hipError_t launch2_col(int op, int grid, const Col2Args& a, hipStream_t s);
template <int H>
hipError_t launch2_row(int mode, int grid, const Row2Args& a, hipStream_t s);

// direct (FFT-free) A x (transpose = 0) or A^T r (transpose = 1), d in
// {2, 4, 8, 16} (inst_direct.hip)
hipError_t launch_direct(int transpose, int d, const float* c, const float* in, float* out, long long n,
                         hipStream_t s);

}  // namespace cs
