// zmc_rtc.hpp -- run-time compiled user integrands (see zmc_rtc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "zmc_device.hpp"

namespace zmc {

constexpr int kUserBase = 100;          // ids of user integrands start here
constexpr int kMaxUserIntegrands = 64;

// Register a body; compiles it once to check it.  ZMC_EINVAL with the
// compiler log in the thread's error text when it does not compile.
int rtc_register(const char* body, int n_params, int* id);
// n_params of a registered user integrand, -1 if unknown.
int rtc_n_params(int id);
// Launch the (id, dim, eval) sampling kernel (compiled on first use) over
// the a.total_units units from a.unit0 on, with a persistent grid.
int rtc_launch(int id, int dim, int eval, hipStream_t st, const SampleArgs& a);

} // namespace zmc
