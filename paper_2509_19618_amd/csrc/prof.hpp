// prof.hpp -- optional per-kernel-class timing with HIP events, recorded on
// the stream each kernel is launched on.  Off by default; when on, every
// instrumented launch is bracketed by two events from a reusable pool and
// the elapsed times are folded in when the caller collects (after it has
// synchronised the stream).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mxp {
namespace prof {

enum Cls : int { GEMM = 0, TRSM = 1, DIAG = 2, PREC = 3, REGEN = 4, GMRES = 5, GEMM64 = 6, NCLS = 7 };

bool enabled();
// begin() records a start event on s and returns it (nullptr when timing of
// class c is off); end() records the matching stop event on the same stream.
hipEvent_t begin(Cls c, hipStream_t s);
void end(hipEvent_t start, Cls c, hipStream_t s, double flops, double bytes);

}  // namespace prof
}  // namespace mxp
