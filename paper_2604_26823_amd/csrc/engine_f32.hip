// FP32 instantiation of the hot-path engine.
#include "engine_impl.h"

namespace ic {
template <>
size_t workspace_bytes_t<float>(const ic_problem& p) {
  Engine<float> e(p, nullptr, 0, nullptr);
  return e.needed();
}
template <>
EngineBase* make_engine_t<float>(const ic_problem& p, void* ws, size_t ws_bytes,
                                 hipStream_t stream) {
  return new Engine<float>(p, static_cast<char*>(ws), ws_bytes, stream);
}
}  // namespace ic
