// C entry points of the batched compression (include/rsvd.h) and the HIP
// graph wrapper used to replay it.
#include <new>

#include "../../include/rsvd.h"
#include "internal.hpp"

using namespace rsvd;

namespace {

inline size_t rup(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct BatchedLayout {
  size_t order, queue, scratch, total;
};

BatchedLayout batched_layout(int nblk, int nwg) {
  BatchedLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off = rup(off + b, 256); return o; };
  L.order = take((size_t)nblk * sizeof(int));
  L.queue = take(256);
  L.scratch = take((size_t)nwg * batched_scratch_doubles_per_wg() * sizeof(double));
  L.total = off;
  return L;
}

int default_wg() {
  int dev = 0, cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      cu = prop.multiProcessorCount;
  }
  return 2 * cu;
}

}  // namespace

struct rsvd_graph_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

rsvd_status rsvd_batched_workspace_size(int32_t nblk, int32_t n_workgroups, size_t* h_bytes) {
  if (!h_bytes || nblk < 1 || n_workgroups < 0 || n_workgroups > 65536) return RSVD_E_ARG;
  int nwg = n_workgroups ? n_workgroups : default_wg();
  *h_bytes = batched_layout(nblk, nwg).total;
  return RSVD_OK;
}

rsvd_status rsvd_batched(int32_t nblk, const int32_t* d_m, const int32_t* d_n, const float* const* d_A,
                         const int32_t* d_lda, double eps, int32_t rank_cap, uint64_t seed, float* d_U, double* d_S,
                         float* d_V, const int64_t* d_offU, const int64_t* d_offV, int32_t* d_rank,
                         int32_t* d_status, int32_t n_workgroups, void* d_ws, size_t ws_bytes, void* stream) {
  if (nblk < 1 || !d_m || !d_n || !d_A || !d_lda || !d_U || !d_S || !d_V || !d_offU || !d_offV || !d_rank ||
      !d_status)
    return RSVD_E_ARG;
  if (!(eps > 0.0) || !(eps < 1.0) || rank_cap < 16 || rank_cap > batched_max_rank() || n_workgroups < 0 ||
      n_workgroups > 65536)
    return RSVD_E_ARG;
  int nwg = n_workgroups ? n_workgroups : default_wg();
  BatchedLayout L = batched_layout(nblk, nwg);
  if (!d_ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return RSVD_E_WORKSPACE;
  char* ws = reinterpret_cast<char*>(d_ws);
  hipError_t e = launch_batched(nblk, d_m, d_n, d_A, d_lda, eps, rank_cap, seed, d_U, d_S, d_V, d_offU, d_offV,
                                d_rank, d_status, reinterpret_cast<int*>(ws + L.order),
                                reinterpret_cast<int*>(ws + L.queue), reinterpret_cast<double*>(ws + L.scratch), nwg,
                                reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? RSVD_OK : RSVD_E_HIP;
}

rsvd_status rsvd_batched_graph_create(int32_t nblk, const int32_t* d_m, const int32_t* d_n,
                                      const float* const* d_A, const int32_t* d_lda, double eps, int32_t rank_cap,
                                      uint64_t seed, float* d_U, double* d_S, float* d_V, const int64_t* d_offU,
                                      const int64_t* d_offV, int32_t* d_rank, int32_t* d_status,
                                      int32_t n_workgroups, void* d_ws, size_t ws_bytes, void* stream,
                                      rsvd_graph_t* h_out) {
  if (!h_out) return RSVD_E_ARG;
  *h_out = nullptr;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (st == nullptr) return RSVD_E_ARG;   // the legacy default stream cannot be captured
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return RSVD_E_HIP;
  rsvd_status s = rsvd_batched(nblk, d_m, d_n, d_A, d_lda, eps, rank_cap, seed, d_U, d_S, d_V, d_offU, d_offV,
                               d_rank, d_status, n_workgroups, d_ws, ws_bytes, stream);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(st, &graph);
  if (s != RSVD_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess || !graph) return RSVD_E_HIP;
  rsvd_graph_s* g = new (std::nothrow) rsvd_graph_s();
  if (!g) { (void)hipGraphDestroy(graph); return RSVD_E_HIP; }
  g->graph = graph;
  if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    delete g;
    return RSVD_E_HIP;
  }
  *h_out = g;
  return RSVD_OK;
}

rsvd_status rsvd_graph_launch(rsvd_graph_t g, void* stream) {
  if (!g) return RSVD_E_ARG;
  return hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? RSVD_OK : RSVD_E_HIP;
}

void rsvd_graph_destroy(rsvd_graph_t g) {
  if (!g) return;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
