// A captured cycle: the launches of one cycle recorded once into a HIP graph
// and replayed once per cycle.
#pragma once
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "h2_impl.h"

namespace h2mg {

struct CycleGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  CycleGraph() = default;
  CycleGraph(const CycleGraph&) = delete;
  CycleGraph& operator=(const CycleGraph&) = delete;
  ~CycleGraph() { reset(); }
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};

// Record the launches of body() into g on the handle's private capture
// stream (the caller's stream may be the null stream, which cannot be
// captured), then instantiate it.
template <typename F>
void capture(H2& h, CycleGraph& g, F&& body) {
  auto check = [](hipError_t e, const char* what) {
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
  };
  hipStream_t user = h.stream;
  if (!h.capture_stream) check(hipStreamCreateWithFlags(&h.capture_stream, hipStreamNonBlocking), "stream create");
  h.stream = h.capture_stream;
  check(hipStreamBeginCapture(h.capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  try {
    body();
  } catch (...) {
    hipGraph_t partial = nullptr;
    (void)hipStreamEndCapture(h.capture_stream, &partial);
    if (partial) (void)hipGraphDestroy(partial);
    h.stream = user;
    throw;
  }
  h.stream = user;
  check(hipStreamEndCapture(h.capture_stream, &g.graph), "end capture");
  check(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0), "graph instantiate");
}

}  // namespace h2mg
