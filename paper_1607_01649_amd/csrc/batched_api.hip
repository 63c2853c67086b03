// C entry points of the batched compression (include/rsvd.h) and the HIP
// graph wrapper used to replay it.
#include <algorithm>
#include <new>
#include <vector>

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

// One persistent workgroup per resident slot: compute units x workgroups that fit on one.
int default_wg() {
  int dev = 0, cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      cu = prop.multiProcessorCount;
  }
  return cu * batched_resident_per_cu();
}

bool tiles_valid(const int32_t* t) {
  if (!t) return true;
  for (int c = 0; c < RSVD_BATCHED_CLASSES; ++c)
    if (t[c] < 0 || t[c] >= RSVD_BATCHED_TILE_VARIANTS) return false;
  return true;
}

struct BatchedCall {
  int32_t nblk;
  const int32_t *m, *n;
  const float* const* A;
  const int32_t* lda;
  double eps;
  int32_t rank_cap;
  uint64_t seed;
  float* U;
  double* S;
  float* V;
  const int64_t *offU, *offV;
  int32_t *rank, *status;
  int32_t n_workgroups;
  void* ws;
  size_t ws_bytes;
};

rsvd_status batched_check(const BatchedCall& c) {
  if (c.nblk < 1 || !c.m || !c.n || !c.A || !c.lda || !c.U || !c.S || !c.V || !c.offU || !c.offV || !c.rank ||
      !c.status)
    return RSVD_E_ARG;
  if (!(c.eps > 0.0) || !(c.eps < 1.0) || c.rank_cap < 16 || c.rank_cap > batched_max_rank() ||
      c.n_workgroups < 0 || c.n_workgroups > 65536)
    return RSVD_E_ARG;
  const int nwg = c.n_workgroups ? c.n_workgroups : default_wg();
  if (!c.ws || c.ws_bytes < batched_layout(c.nblk, nwg).total || (reinterpret_cast<uintptr_t>(c.ws) & 255) != 0)
    return RSVD_E_WORKSPACE;
  return RSVD_OK;
}

hipError_t batched_launch(const BatchedCall& c, const int* tiles, int class_mask, hipStream_t st) {
  const int nwg = c.n_workgroups ? c.n_workgroups : default_wg();
  const BatchedLayout L = batched_layout(c.nblk, nwg);
  char* ws = reinterpret_cast<char*>(c.ws);
  return launch_batched(c.nblk, c.m, c.n, c.A, c.lda, c.eps, c.rank_cap, c.seed, c.U, c.S, c.V, c.offU, c.offV,
                        c.rank, c.status, reinterpret_cast<int*>(ws + L.order), reinterpret_cast<int*>(ws + L.queue),
                        reinterpret_cast<double*>(ws + L.scratch), nwg, tiles, class_mask, st);
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
                         int32_t* d_status, int32_t n_workgroups, const int32_t* h_tiles, void* d_ws,
                         size_t ws_bytes, void* stream) {
  const BatchedCall c{nblk, d_m, d_n, d_A, d_lda, eps, rank_cap, seed, d_U, d_S, d_V, d_offU, d_offV,
                      d_rank, d_status, n_workgroups, d_ws, ws_bytes};
  const rsvd_status s = batched_check(c);
  if (s != RSVD_OK) return s;
  if (!tiles_valid(h_tiles)) return RSVD_E_ARG;
  return batched_launch(c, h_tiles, (1 << RSVD_BATCHED_CLASSES) - 1, reinterpret_cast<hipStream_t>(stream)) ==
                 hipSuccess
             ? RSVD_OK
             : RSVD_E_HIP;
}

rsvd_status rsvd_batched_autotune(int32_t nblk, const int32_t* d_m, const int32_t* d_n, const float* const* d_A,
                                  const int32_t* d_lda, double eps, int32_t rank_cap, uint64_t seed, float* d_U,
                                  double* d_S, float* d_V, const int64_t* d_offU, const int64_t* d_offV,
                                  int32_t* d_rank, int32_t* d_status, int32_t n_workgroups, void* d_ws,
                                  size_t ws_bytes, void* stream, int32_t* h_tiles_out, float* h_ms_out) {
  if (!h_tiles_out) return RSVD_E_ARG;
  const BatchedCall c{nblk, d_m, d_n, d_A, d_lda, eps, rank_cap, seed, d_U, d_S, d_V, d_offU, d_offV,
                      d_rank, d_status, n_workgroups, d_ws, ws_bytes};
  rsvd_status s = batched_check(c);
  if (s != RSVD_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  constexpr int NC = RSVD_BATCHED_CLASSES, NV = RSVD_BATCHED_TILE_VARIANTS;
  const int def = batched_default_variant();
  // blocks per size class (the same classes the kernel uses: max(m, n) in 128-wide bins)
  std::vector<int32_t> hm(nblk), hn(nblk);
  if (hipMemcpyAsync(hm.data(), d_m, sizeof(int32_t) * nblk, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(hn.data(), d_n, sizeof(int32_t) * nblk, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return RSVD_E_HIP;
  int count[NC] = {0};
  for (int b = 0; b < nblk; ++b) {
    const int mx = std::max(hm[b], hn[b]);
    if (mx >= 1 && mx <= batched_max_dim()) ++count[(mx - 1) >> 7];
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return RSVD_E_HIP;
  }
  constexpr int kReps = 2;
  int tiles[NC];
  for (int k = 0; k < NC; ++k) tiles[k] = def;
  s = RSVD_OK;
  for (int cls = 0; cls < NC && s == RSVD_OK; ++cls) {
    float best = 0.f;
    int bestv = def;
    for (int v = 0; v < NV && s == RSVD_OK; ++v) {
      float ms = 0.f;
      if (count[cls] > 0) {
        int trial[NC];
        for (int k = 0; k < NC; ++k) trial[k] = def;
        trial[cls] = v;
        bool ok = batched_launch(c, trial, 1 << cls, st) == hipSuccess;   // warm-up
        ok = ok && hipEventRecord(e0, st) == hipSuccess;
        for (int r = 0; r < kReps && ok; ++r) ok = batched_launch(c, trial, 1 << cls, st) == hipSuccess;
        ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (!ok) { s = RSVD_E_HIP; break; }
        ms /= kReps;
        if (v == 0 || ms < best) { best = ms; bestv = v; }
      }
      if (h_ms_out) h_ms_out[cls * NV + v] = ms;
    }
    tiles[cls] = bestv;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != RSVD_OK) return s;
  for (int k = 0; k < NC; ++k) h_tiles_out[k] = tiles[k];
  return RSVD_OK;
}

rsvd_status rsvd_batched_graph_create(int32_t nblk, const int32_t* d_m, const int32_t* d_n,
                                      const float* const* d_A, const int32_t* d_lda, double eps, int32_t rank_cap,
                                      uint64_t seed, float* d_U, double* d_S, float* d_V, const int64_t* d_offU,
                                      const int64_t* d_offV, int32_t* d_rank, int32_t* d_status,
                                      int32_t n_workgroups, const int32_t* h_tiles, void* d_ws, size_t ws_bytes,
                                      void* stream, rsvd_graph_t* h_out) {
  if (!h_out) return RSVD_E_ARG;
  *h_out = nullptr;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (st == nullptr) return RSVD_E_ARG;   // the legacy default stream cannot be captured
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return RSVD_E_HIP;
  rsvd_status s = rsvd_batched(nblk, d_m, d_n, d_A, d_lda, eps, rank_cap, seed, d_U, d_S, d_V, d_offU, d_offV,
                               d_rank, d_status, n_workgroups, h_tiles, d_ws, ws_bytes, stream);
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
