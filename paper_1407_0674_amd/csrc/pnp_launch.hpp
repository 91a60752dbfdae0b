// The launch table of the evaluation's passes for one (precision, grid
// size, launch variant): host functions that launch each pass kernel over a
// device table of per-instance arguments.  The tables of each (precision,
// size, FFT schedule) are built in their own translation unit (pnp_ops.hip
// compiled once per triple), so they compile in parallel; the ABI's
// translation unit only declares ops_inst.
#pragma once
#include <hip/hip_runtime.h>

#include "pnp_kernels.hpp"

namespace pnp {

struct Ops {
  void (*tables)(const TableArgs*, int, int, int, hipStream_t);
  void (*zfwd)(const EvalArgs*, int, hipStream_t);
  void (*ystep)(const EvalArgs*, int, int, int, bool, int, hipStream_t);  // count, sel, nf, fwd, part
  void (*xfwd)(const EvalArgs*, int, int, hipStream_t);                   // count, part
  void (*zderiv)(const EvalArgs*, int, bool, int, hipStream_t);
  void (*xback)(const EvalArgs*, int, int, bool, int, hipStream_t);  // count, smax, large, part
  int zderiv_tiles;  // workgroups of the derivative pass per instance
  void (*zinv)(const EvalArgs*, int, int, hipStream_t);
  void (*xplain)(const EvalArgs*, int, int, bool, hipStream_t);
  void (*xport)(const EvalArgs*, int, double*, int, hipStream_t);
  uint32_t sched_alt;  // passes (bit p: pass p) whose secondary FFT schedule differs from the primary
};

// Grids up to kNarrowMax also have the narrow tile shape (V bit 0); larger
// ones already launch thousands of workgroups per pass.  Every size has both
// FFT schedules (V bit 1).
constexpr int kNarrowMax = 128;

// the launch table of (T, N, V); defined by the translation unit of
// (T, N, schedule)
template <typename T, int N, int V> const Ops* ops_inst();

}  // namespace pnp
