// Checked kernel launch, used by the launcher sections of the kernel files.
#pragma once

#include "dtw_internal.h"

namespace dtw {

// Launch `fn` on `st` after check_launch has accepted the configuration; the
// arguments are converted to the kernel's parameter types.
template <typename... P, typename... A>
hipError_t launch_checked(void (*fn)(P...), int grid, int threads, size_t dyn_lds, hipStream_t st, A&&... args) {
  const hipError_t e = check_launch(reinterpret_cast<const void*>(fn), grid, threads, dyn_lds);
  if (e != hipSuccess) return e;
  fn<<<grid, threads, dyn_lds, st>>>(static_cast<P>(args)...);
  return hipGetLastError();
}

}  // namespace dtw
