// One path for the kernel launches of the aggregator forward: straight onto a
// stream, or, while a Recording is active on the calling thread, into that
// recording (the graph mode of the aggregate entry points replays recordings
// as HIP graphs).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <tuple>
#include <utility>
#include <vector>

namespace vggtx {

// One recorded launch: the kernel, its shape and its argument bytes (each
// argument at an offset aligned for its type, padding zeroed).
struct LaunchRecord {
  const void* func = nullptr;
  dim3 grid, block;
  unsigned shm = 0;
  std::vector<uint8_t> args;
  std::vector<uint32_t> offs;
};

struct Recording {
  std::vector<LaunchRecord> launches;
};

// The recording of the calling thread, or null (launch immediately).
Recording*& active_recording();

namespace detail {
template <typename Tuple, size_t... I>
hipError_t launch_now(const void* f, dim3 g, dim3 b, unsigned shm, hipStream_t s, Tuple& t,
                      std::index_sequence<I...>) {
  void* argv[] = {(void*)&std::get<I>(t)..., nullptr};
  return hipLaunchKernel(f, g, b, argv, shm, s);
}

template <typename Tuple, size_t... I>
void record(const void* f, dim3 g, dim3 b, unsigned shm, Tuple& t, std::index_sequence<I...>) {
  LaunchRecord r;
  r.func = f;
  r.grid = g;
  r.block = b;
  r.shm = shm;
  size_t off = 0;
  auto put = [&](const auto& v) {
    const size_t al = alignof(std::decay_t<decltype(v)>);
    off = (off + al - 1) / al * al;
    r.offs.push_back((uint32_t)off);
    if (r.args.size() < off + sizeof(v)) r.args.resize(off + sizeof(v), 0);
    memcpy(r.args.data() + off, &v, sizeof(v));
    off += sizeof(v);
  };
  (put(std::get<I>(t)), ...);
  active_recording()->launches.push_back(std::move(r));
}
}  // namespace detail

// Launch `kernel` with the arguments converted to its parameter types.
template <typename... P, typename... A>
hipError_t launch(void (*kernel)(P...), dim3 grid, dim3 block, unsigned shm, hipStream_t s, A&&... a) {
  static_assert(sizeof...(P) == sizeof...(A), "argument count");
  std::tuple<P...> t(static_cast<P>(std::forward<A>(a))...);
  if (active_recording()) {
    detail::record((const void*)kernel, grid, block, shm, t, std::index_sequence_for<P...>{});
    return hipSuccess;
  }
  return detail::launch_now((const void*)kernel, grid, block, shm, s, t, std::index_sequence_for<P...>{});
}

}  // namespace vggtx
