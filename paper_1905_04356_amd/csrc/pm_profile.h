// pm_profile.h -- optional per-kernel device timing with HIP events, and the
// launch helper every kernel of the library goes through.
#pragma once
#include <hip/hip_runtime.h>

#include <tuple>
#include <type_traits>
#include <utility>

namespace pm {

enum KernelKind {
  K_NTT_FWD = 0, K_POINTWISE = 1, K_NTT_INV = 2, K_CRT = 3, K_BATCHED = 4,
  K_VDM_EVAL = 5, K_VDM_INTERP = 6, K_GEO = 7
};

bool profiling();

// A timing scope.  By default launches made through launch() inside it are
// timed as `kind`, each by events that its own dispatch fills, which puts no
// extra packets on the stream.  With scope_events the whole scope is timed
// by an event pair instead: for graph replays, whose kernels do not pass
// through launch().  Nothing is timed inside a stream capture.
class KernelTimer {
 public:
  KernelTimer(int kind, hipStream_t s, bool scope_events = false);
  ~KernelTimer();
  KernelTimer(const KernelTimer&) = delete;
  KernelTimer& operator=(const KernelTimer&) = delete;

 private:
  int kind_;
  int prev_kind_;
  hipStream_t s_;
  hipEvent_t a_{}, b_{};
  bool armed_ = false;
};

// Launch the kernel at `fn` with argument pointers `args`; returns the
// launch's error, else the last error HIP holds (which it clears).
hipError_t launch_kernel(const void* fn, dim3 grid, dim3 block, void** args, size_t lds,
                         hipStream_t s);

namespace detail {
template <typename Tuple, size_t... I>
void arg_ptrs(Tuple& t, void** p, std::index_sequence<I...>) {
  ((p[I] = (void*)&std::get<I>(t)), ...);
}
}  // namespace detail

// Typed form: converts the arguments to the kernel's parameter types.
template <typename... Params, typename... Args>
hipError_t launch(void (*kernel)(Params...), dim3 grid, dim3 block, size_t lds, hipStream_t s,
                  Args&&... args) {
  static_assert(sizeof...(Params) == sizeof...(Args), "kernel argument count");
  std::tuple<std::decay_t<Params>...> vals{std::forward<Args>(args)...};
  void* ptrs[sizeof...(Params) > 0 ? sizeof...(Params) : 1];
  detail::arg_ptrs(vals, ptrs, std::index_sequence_for<Params...>{});
  return launch_kernel((const void*)kernel, grid, block, ptrs, lds, s);
}

}  // namespace pm
